"""Adaptive Dormand-Prince 5(4) stepping on the GPU against the oracle.

Two instances (Schwarzschild and spin 0.5) advance one attempt at a time with
their own steps; the first is perturbed and starts with an overlong step, so
it is rejected before it is accepted.  Every attempt is checked from the same
inputs on both sides (the GPU's state, steps and rejection flags before it):
identical accept decisions and a state equal to the oracle's to 1e-12 of its
scale.  The error norm and the next step are compared to 1e-6 relative: the
norm measures the difference of the fifth- and fourth-order solutions, which
near the tolerance is about 1e-5 of the step's change dt |L(u)|, so the
1e-12 relative parity of the stage derivatives leaves it about 1e-7 relative
(the next step follows it through err^-1/5).
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain, dp5  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def _setup(shells, holes, filt, pert_amp=1e-2):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = len(holes)
    wl = configs.Workload("dp5", shells, holes, [(1.0, -1.0, 1.0)] * n, [0.01] * n, filt, 1, None)
    d = domain.Domain([domain.Shell(*s) for s in shells], filter_params=filt)
    u0, ubg, H, dH = wl.initial_data(d.xyz(), d.offsets)
    owner = d.instance_of_value()
    u0 = u0 + np.where(owner == 0, d.to_layout(inputs.smooth_random_field(d.xyz(), pert_amp, 3, 3, 2.0)), 0.0)
    s = ghmi.GHSolver(shells, n, filt)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    return wl, d, s, u0, ubg, H, dH


SHELLS = [(0, 7, 5, 1.8, 3.0), (0, 7, 5, 3.0, 4.5), (1, 7, 3, 1.7, 3.2)]
HOLES = [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0, 0, 1))]


def _run(wl, d, s, u0, ubg, H, dH, dt0, atol, rtol, n):
    u = dev(u0)
    t = torch.zeros(wl.n_inst, dtype=torch.float64, device="cuda:0")
    dt = dev(np.array(dt0, dtype=float))
    rej = torch.zeros(wl.n_inst, dtype=torch.int32, device="cuda:0")
    na = torch.zeros(wl.n_inst, dtype=torch.int32, device="cuda:0")
    err = torch.zeros(wl.n_inst, dtype=torch.float64, device="cuda:0")
    n_rej = 0
    for a in range(n):
        u_in, dt_in, rej_in = u.cpu().numpy(), dt.cpu().numpy(), rej.cpu().numpy().astype(bool)
        t_in, na_in = t.cpu().numpy(), na.cpu().numpy()
        s.step_dp5(u, 1, atol, rtol, t, dt, rejected=rej, n_accepted=na, err=err)
        acc_g = (na.cpu().numpy() - na_in) > 0
        uo, acc_o, dt_o, err_o = d.dp5_attempt(u_in, H, dH, ubg, wl.gamma, dt_in, atol, rtol, rej_in)
        n_rej += int((~acc_o).sum())
        assert np.array_equal(acc_g, acc_o), (a, acc_g, acc_o, err.cpu().numpy(), err_o)
        assert np.array_equal(rej.cpu().numpy().astype(bool), ~acc_o)
        assert np.allclose(err.cpu().numpy(), err_o, rtol=1e-6, atol=0), (a, err.cpu().numpy(), err_o)
        assert np.allclose(dt.cpu().numpy(), dt_o, rtol=1e-6, atol=0), (a, dt.cpu().numpy(), dt_o)
        assert np.array_equal(t.cpu().numpy(), t_in + np.where(acc_o, dt_in, 0.0))
        diff = np.max(np.abs(u.cpu().numpy() - uo))
        assert diff <= 1e-12 * np.max(np.abs(uo)), (a, diff)
    return n_rej, t.cpu().numpy(), dt.cpu().numpy()


def test_dp5_attempts_match_oracle_with_rejections():
    wl, d, s, u0, ubg, H, dH = _setup(SHELLS, HOLES, None)
    n_rej, t, dt = _run(wl, d, s, u0, ubg, H, dH, [0.3, 0.02], 1e-8, 1e-8, 8)
    print(f"  8 attempts: {n_rej} rejections, t = {t}, dt = {dt}", flush=True)
    assert n_rej >= 1 and np.all(t > 0)


def test_dp5_with_filter_matches_oracle():
    rs = configs.geometric_radii(1.8, 6.0, 2)
    shells = [(0, 9, 7, rs[0], rs[1]), (0, 9, 7, rs[1], rs[2])]
    wl, d, s, u0, ubg, H, dH = _setup(shells, [(1.0, 0.3, (0.2, 0.1, 1.0))], configs.FILTER_DEFAULT, 1e-3)
    n_rej, t, dt = _run(wl, d, s, u0, ubg, H, dH, [0.05], 1e-9, 1e-9, 6)
    print(f"  6 filtered attempts: {n_rej} rejections, t = {t}", flush=True)
    assert t[0] > 0


def test_one_call_of_n_attempts_equals_n_calls():
    """The first-same-as-last reuse inside one call gives bitwise the state of
    separate calls (which evaluate the first stage anew) that pass the
    rejection flags on."""
    wl, d, s, u0, ubg, H, dH = _setup(SHELLS, HOLES, None, 1e-4)
    outs = []
    for calls in ((4,), (1, 1, 1, 1)):
        u = dev(u0)
        t = torch.zeros(2, dtype=torch.float64, device="cuda:0")
        dt = dev(np.array([0.002, 0.002]))
        na = torch.zeros(2, dtype=torch.int32, device="cuda:0")
        rej = torch.zeros(2, dtype=torch.int32, device="cuda:0")
        for n in calls:
            s.step_dp5(u, n, 1e-6, 1e-6, t, dt, rejected=rej, n_accepted=na)
        assert na.cpu().tolist() == [4, 4]
        outs.append((u, t, dt))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_dp5_argument_errors():
    wl, d, s, u0, ubg, H, dH = _setup(SHELLS, HOLES, None)
    u = dev(u0)
    t = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    dt = dev(np.array([0.01, 0.01]))
    for bad in ((-1, 1e-8, 1e-8), (1, 0.0, 0.0), (1, -1e-8, 1e-8), (1, float("nan"), 1e-8)):
        with pytest.raises(ghmi.GHError) as ei:
            s.step_dp5(u, bad[0], bad[1], bad[2], t, dt)
        assert ei.value.code == -1
    assert dp5.MINSCALE == 0.2

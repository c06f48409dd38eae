"""The workloads at their stated lengths, and the two-level checkpoint
schedule of the reverse pass on the GPU.

* The 8-shell pulse workload for its 1000 RK3 steps and the 20-shell L = 31
  domain for its 2000 (unfiltered): the state stays finite, and the
  constraint norm stays bounded (the damped system keeps it from growing).
  The 20-shell run answers the question whether unfiltered evolutions drift
  through the half of the angular grid values the Y_lm derivatives do not
  see: if they did, the norm would grow and a projection after every step
  would be needed.
* A two-level schedule (inner checkpoints inside each outer segment) gives
  bitwise the gradient of the one-level schedule: the recomputed states are
  the same deterministic steps.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_1804_09101_amd import autograd as gha  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _upload(wl):
    xyz = ghmi.grid_coords(wl.shells)
    offs = np.concatenate([[0], np.cumsum([s[1] * 2 * (s[2] + 1) ** 2 for s in wl.shells])])
    u0, ubg, H, dH = wl.initial_data(xyz, offs, device="cuda:0")
    s = ghmi.GHSolver(wl.shells, wl.n_inst, wl.filter_params)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    return s, dev(u0)


def _norm(s, u):
    return float(s.constraints(u, want_C=False)[1].cpu()[0])


def test_pulse_8shell_1000_steps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = configs.pulse_8shell()
    print(f"\n[case] pulse_8shell, {wl.n_steps} RK3 steps", flush=True)
    s, u0 = _upload(wl)
    u = u0.clone()
    n0 = _norm(s, u)
    norms = []
    for _ in range(4):
        s.step(u, wl.n_steps // 4)
        norms.append(_norm(s, u))
        print(f"  constraint norm {norms[-1]:.3e} (start {n0:.3e})", flush=True)
    assert bool(torch.isfinite(u).all())
    change = float((u - u0).abs().max())
    print(f"  max change {change:.3e}", flush=True)
    assert max(norms) < 2.0 * n0 and change < 1e-2
    s.close()


def test_large_20shell_2000_steps_unfiltered():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = configs.large_20shell()
    print(f"\n[case] large_20shell, {wl.n_steps} RK3 steps, no filter", flush=True)
    s, u0 = _upload(wl)
    s.set_angular(2)               # the faster form of the same operators
    u = u0.clone()
    n0 = _norm(s, u)
    norms = []
    for _ in range(8):
        s.step(u, wl.n_steps // 8)
        norms.append(_norm(s, u))
        print(f"  constraint norm {norms[-1]:.3e} (start {n0:.3e})", flush=True)
    assert bool(torch.isfinite(u).all())
    change = float((u - u0).abs().max())
    print(f"  max change {change:.3e}", flush=True)
    assert max(norms) < 2.0 * n0 and change < 1e-3
    s.close()


def test_two_level_schedule_gives_the_one_level_gradient():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rs = configs.geometric_radii(1.8, 6.0, 2)
    shells = [(0, 9, 5, rs[0], rs[1]), (0, 9, 5, rs[1], rs[2])]
    wl = configs.Workload("ckpt", shells, [(1.0, 0.3, (0, 0, 1))], [(0.9, -0.5, 1.2)], [0.006],
                          configs.FILTER_DEFAULT, 1, None)
    print("\n[case] two-level checkpoints: 24 steps, k = 8 against k1 = 12, k2 = 3", flush=True)
    s, u0 = _upload(wl)
    xyz = ghmi.grid_coords(shells)
    offs = np.concatenate([[0], np.cumsum([sh[1] * 2 * (sh[2] + 1) ** 2 for sh in shells])])
    u0 = u0 + dev(configs.to_layout(inputs.smooth_random_field(xyz, 1e-2, 3, 3, 2.0), shells, offs))
    grads = []
    for k1, k2 in ((8, None), (12, 3), (24, 5)):
        gamma = torch.tensor(wl.gamma, dtype=torch.float64, requires_grad=True)
        ua = u0.clone().requires_grad_(True)
        un = gha.evolve(ua, gamma, s, wl.dt, 24, checkpoint_every=k1, save_derivatives=False, inner_every=k2)
        gha.constraint_norm(un, s).sum().backward()
        grads.append((ua.grad.clone(), gamma.grad.clone()))
    for gu, gg in grads[1:]:
        assert torch.equal(gu, grads[0][0]) and torch.equal(gg, grads[0][1])
    assert float(grads[0][0].abs().max()) > 0
    s.close()

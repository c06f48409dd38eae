"""The SSP-RK3 stages of a step against gh_rhs on the stage states.

In a step the pointwise kernel writes the new state of every point off the
treated faces itself, and a face kernel applies the boundary treatment to the
interface and outer faces and finishes them; gh_rhs instead writes d_t u
everywhere and treats the faces with its own boundary kernel.  So each stage
that gh_step_stages stores must equal c0 u0 + c1 (us + dt gh_rhs(us)) to
rounding: stage 1 with (c0, c1) = (0, 1), stage 2 (3/4, 1/4), stage 3 (1/3,
2/3), for every combination of the outer boundary (Dirichlet or
constraint-preserving) and of the interface projection (frozen or from the
state), on two instances with interfaces and per-instance time steps.  A wrong
face set or a missed stage term moves the state by O(dt |L|), about 1e-3 of
its size here; the bar is 1e-13 of the state.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu

SHELLS = [(0, 9, 7, 1.8, 3.0), (0, 9, 7, 3.0, 4.6), (0, 8, 7, 4.6, 6.0),
          (1, 7, 5, 1.5, 2.9), (1, 9, 5, 2.9, 5.0)]
HOLES = [(1.0, 0.0, (0.0, 0.0, 1.0)), (0.9, 0.5, (0.3, -0.2, 0.9))]
GAMMA = [(1.0, 0.5, 1.0), (0.7, -1.0, 1.3)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def test_step_stages_equal_rhs_stage_updates():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dt = [configs.COURANT * min(configs.min_radial_spacing(s[1], s[3], s[4]) for s in SHELLS if s[0] == i)
          for i in range(2)]
    wl = configs.Workload("stage_split", SHELLS, HOLES, GAMMA, dt, None, 1, None)
    xyz = ghmi.grid_coords(SHELLS)
    offs = np.concatenate([[0], np.cumsum([s[1] * 2 * (s[2] + 1) ** 2 for s in SHELLS])])
    u0, ubg, H, dH = wl.initial_data(xyz, offs)
    u0 = u0 + configs.to_layout(inputs.smooth_random_field(xyz, 1e-2, 5, 3, 2.0), SHELLS, offs)
    # the time step of each field element: its shell's instance's
    dtf = dev(np.concatenate([np.full(50 * (offs[k + 1] - offs[k]), dt[sh[0]]) for k, sh in enumerate(SHELLS)]))
    u = dev(u0)
    scale = float(u.abs().max())
    finals = {}
    for outer_mode in (0, 1):
        for iface_mode in (0, 1):
            print(f"\n[case] stage split: outer_mode {outer_mode}, interface mode {iface_mode}", flush=True)
            s = ghmi.GHSolver(SHELLS, 2, None)
            s.set_background(dev(H), dev(dH), dev(ubg))
            s.set_params(wl.gamma, wl.dt)
            s.set_outer_bc(outer_mode)
            s.set_interface(iface_mode)
            un = u.clone()
            u1, u2 = torch.empty_like(u), torch.empty_like(u)
            s.step_stages(un, u1, u2)
            stages = ((0.0, 1.0, u, u1), (0.75, 0.25, u1, u2), (1.0 / 3.0, 2.0 / 3.0, u2, un))
            for k, (c0, c1, us, got) in enumerate(stages):
                ref = c1 * (us + dtf * s.rhs(us))
                if c0:
                    ref = ref + c0 * u
                err = float((got - ref).abs().max()) / scale
                moved = float((got - us).abs().max()) / scale
                print(f"  stage {k + 1}: |step stage - rhs stage| {err:.2e} of the state (the stage moves it by "
                      f"{moved:.1e})", flush=True)
                assert err < 1e-13 and moved > 1e-6
            finals[(outer_mode, iface_mode)] = un
            s.close()
    # both switches change the step (so both face paths ran)
    d_outer = float((finals[(1, 0)] - finals[(0, 0)]).abs().max()) / scale
    d_iface = float((finals[(0, 1)] - finals[(0, 0)]).abs().max()) / scale
    print(f"  step difference: outer mode {d_outer:.2e}, interface mode {d_iface:.2e} of the state", flush=True)
    assert d_outer > 1e-12 and d_iface > 1e-14

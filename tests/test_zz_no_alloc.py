"""gh_constraints_static (partial sums in a file-scope device array, no
allocation in the call) against gh_constraints on the same inputs, through the
C interface: the constraints and the norm must be bitwise equal.  Two calls in
a row, the second on a smaller domain (another context on the same GPU, so
the shared array holds the first call's partial sums when it starts)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _case(shells, holes, seed):
    wl = configs.Workload("static", shells, holes, [configs.GAMMA_DEFAULT] * len(holes), [0.005] * len(holes),
                          None, 1, None)
    d = domain.Domain([domain.Shell(*s) for s in shells])
    xyz = d.xyz()
    u0, ubg, H, dH = wl.initial_data(xyz, d.offsets)
    u0 = u0 + d.to_layout(inputs.smooth_random_field(xyz, 1e-2, seed, 3, 2.0))
    s = ghmi.GHSolver(shells, len(holes))
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    return s, dev(u0)


def test_static_scratch_constraints_match_the_allocating_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    big = [(0, 9, 7, 1.8, 3.0), (0, 11, 7, 3.0, 5.0), (1, 7, 5, 1.3, 2.5), (1, 9, 5, 2.5, 4.0)]
    small = [(0, 5, 3, 1.7, 3.0)]
    cases = [(big, [(1.0, 0.3, (0.2, 0.3, 0.9)), (0.8, 0.6, (1.0, 0.0, 0.2))], 1),
             (small, [(1.0, 0.5, (0.0, 0.0, 1.0))], 2)]
    for shells, holes, seed in cases:
        print(f"\n[case] gh_constraints_static, {len(shells)} shells", flush=True)
        s, u = _case(shells, holes, seed)
        C_ref, n_ref = s.constraints(u)
        C = torch.full_like(C_ref, np.nan)
        norm = torch.full_like(n_ref, np.nan)
        torch.cuda.synchronize()
        s.constraints_static(u, C, norm)
        torch.cuda.synchronize()
        print(f"  norm {norm.cpu().numpy()} vs {n_ref.cpu().numpy()}", flush=True)
        assert torch.equal(C, C_ref) and torch.equal(norm, n_ref)
        # the norm alone (no per-point array)
        norm2 = torch.full_like(n_ref, np.nan)
        s.constraints_static(u, None, norm2)
        torch.cuda.synchronize()
        assert torch.equal(norm2, n_ref)
        s.close()

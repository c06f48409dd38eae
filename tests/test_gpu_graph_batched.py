"""Graph replay of whole RK3 steps, and batched instances vs one context per
instance.

* Graph mode replays a captured step; every replay is compared with the eager
  path, with eager torch work and synchronisations between replays.
* A batch of heterogeneous instances in one context (one grouped launch per
  kernel kind) must give exactly the results of one context per instance when
  both run one launch of the same GEMM variant: each output element is then
  accumulated in the same order whatever the tile shape.  With the tuner's
  plans (which may add a tail launch over K chunks, reordering the K sums of
  the last rows) they agree to 1e-13 of the state.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _prepare(wl, pert=1e-3, seed=2):
    d = domain.Domain([domain.Shell(*s) for s in wl.shells], filter_params=wl.filter_params)
    xyz = d.xyz()
    u0, ubg, H, dH = wl.initial_data(xyz, d.offsets)
    u0 = u0 + d.to_layout(inputs.smooth_random_field(xyz, pert, seed, 3, 2.0))
    return d, u0, ubg, H, dH


def _solver(wl, ubg, H, dH):
    s = ghmi.GHSolver(wl.shells, wl.n_inst, wl.filter_params)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    return s


def test_graph_replays_match_eager_steps():
    _need_gpu()
    rs = configs.geometric_radii(1.8, 12.0, 3)
    shells = [(0, 9, 7, rs[i], rs[i + 1]) for i in range(3)]
    wl = configs.Workload("graph", shells, [(1.0, 0.3, (0.2, 0.3, 0.4))], [configs.GAMMA_DEFAULT], [0.004],
                          configs.FILTER_DEFAULT, 1, None)
    d, u0, ubg, H, dH = _prepare(wl)
    eager = _solver(wl, ubg, H, dH)
    graph = _solver(wl, ubg, H, dH)
    graph.set_graph(True)
    ue, ug = dev(u0), dev(u0)
    for chunk in (1, 3, 2, 5):
        eager.step(ue, chunk)
        graph.step(ug, chunk)
        junk = (ug * 2.0).sum() + torch.ones(1000, dtype=torch.float64, device="cuda:0").sum()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert torch.equal(ue, ug), f"graph replay differs after a chunk of {chunk} steps"
    # a new state pointer is captured anew
    ug2 = dev(u0)
    graph.step(ug2, 11)
    torch.cuda.synchronize()
    assert torch.equal(ue, ug2)
    print("  11 steps: graph replays bitwise equal to eager", flush=True)


def test_batched_instances_equal_one_context_per_instance():
    _need_gpu()
    wl = configs.batched_64(seed=3, n_inst=6)
    d, u0, ubg, H, dH = _prepare(wl, pert=1e-4)
    batched = _solver(wl, ubg, H, dH)
    ut = dev(u0)
    batched.step(ut, 3)
    tuned = ut.cpu().numpy()
    pins = [(0, batched.query(6), batched.query(4))]
    if wl.filter_params is not None:
        pins.append((1, batched.query(7), batched.query(5)))
    for p in pins:
        batched.set_gemm_variant(*p)
    ub = dev(u0)
    rhs_b = batched.rhs(ub).cpu().numpy()
    batched.step(ub, 3)
    got = ub.cpu().numpy()
    assert np.max(np.abs(tuned - got)) < 1e-13 * np.max(np.abs(got))
    P = d.P
    for inst in range(wl.n_inst):
        ks = [k for k, s in enumerate(wl.shells) if s[0] == inst]
        sh = [(0,) + tuple(wl.shells[k][1:]) for k in ks]
        lo, hi = 50 * d.offsets[ks[0]], 50 * d.offsets[ks[-1] + 1]
        lo4, hi4 = 4 * d.offsets[ks[0]], 4 * d.offsets[ks[-1] + 1]
        lo16, hi16 = 16 * d.offsets[ks[0]], 16 * d.offsets[ks[-1] + 1]
        wli = configs.Workload("one", sh, [wl.holes[inst]], [wl.gamma[inst]], [wl.dt[inst]], None, 1, None)
        s1 = _solver(wli, ubg[lo:hi], H[lo4:hi4], dH[lo16:hi16])
        for p in pins:
            s1.set_gemm_variant(*p)
        u1 = dev(u0[lo:hi])
        assert np.array_equal(s1.rhs(u1).cpu().numpy(), rhs_b[lo:hi]), inst
        s1.step(u1, 3)
        assert np.array_equal(u1.cpu().numpy(), got[lo:hi]), inst
        s1.close()
    assert P == sum(s[1] * 2 * (s[2] + 1) ** 2 for s in wl.shells)
    print(f"  {wl.n_inst} heterogeneous instances: batched == per-instance, bitwise", flush=True)

"""Every GEMM plan of the library forced into a split plan (gh_set_gemm_plan):
the leading rows in whole rounds of tiles, the remaining rows in smaller tiles
over chunks of K, summed in chunk order.  The autotuner keeps a split only when
it times faster, so these forms are checked here explicitly, with a small
round size so that the test domains' tile counts split.

For each plan the operation that uses it is compared with the oracle at the
usual bars (RHS 1e-12 of the term scale; filters 1e-12 of the state; the
transposes by dot products against the oracle's complex step, 1e-12), and with
the same variant as one launch (the split only reorders the K sums of the
peeled rows: 1e-13)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi, inputs  # noqa: E402

pytestmark = pytest.mark.gpu
H_CS = 1e-30
MIXED = [(0, 9, 7, 1.8, 3.0), (0, 10, 7, 3.0, 5.5), (1, 7, 11, 1.7, 2.9), (1, 6, 11, 2.9, 6.0)]
HOLES = [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0.3, -0.2, 0.9))]
GAMMA = [(0.8, -0.4, 1.2), (1.0, -1.0, 1.0)]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _setup(kind, params):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    wl = configs.Workload("split", MIXED, HOLES, GAMMA, [0.004, 0.004], params, 1, None)
    d = domain.Domain([domain.Shell(*s) for s in MIXED], filter_params=params, filter_kind=kind)
    xyz = d.xyz()
    u0, ubg, H, dH = wl.initial_data(xyz, d.offsets)
    u0 = u0 + d.to_layout(inputs.smooth_random_field(xyz, 1e-2, 5, 3, 2.0))
    s = ghmi.GHSolver(MIXED, 2, params, filter_kind=kind)
    s.set_background(dev(H), dev(dH), dev(ubg))
    s.set_params(wl.gamma, wl.dt)
    return wl, d, s, u0, ubg, H, dH


def _pin_split(s, plan, shape=5):
    """Two K chunks where the tail's K allows (at least 16 per chunk), else one
    (the Fourier GEMMs have K = 2(L+1))."""
    for rnd in (4, 8, 3, 16, 6):
        for chunks in (2, 1):
            try:
                s.set_gemm_plan(plan, shape, 1, 0, chunks, rnd)
                return rnd, chunks
            except ghmi.GHError:
                continue
    raise AssertionError(f"plan {plan}: no round size splits it")


def _term_scale(d, u):
    return max(np.max(np.abs(d.cartesian_derivs(k, b))) for k, b in enumerate(d.split(u, 50)))


def _step_dot(d, s, wl, u0, ubg, H, dH, seed):
    rng = np.random.default_rng(seed)
    lam = rng.standard_normal(u0.shape)
    v = rng.standard_normal(u0.shape)
    jv = d.rk3_step(u0 + 1j * H_CS * v, H, dH, ubg, wl.gamma, wl.dt).imag / H_CS
    ln = s.step_vjp(dev(u0), dev(lam)).cpu().numpy()
    return abs(np.sum(lam * jv) - np.sum(ln * v)) / np.sum(np.abs(lam * jv)), ln


@pytest.mark.parametrize("plan", [0, 1, 2, 3, 4, 5, 6])
def test_split_plans_with_the_exponential_filter(plan):
    wl, d, s, u0, ubg, H, dH = _setup(1, configs.FILTER_DEFAULT)
    print(f"\n[case] forced split of GEMM plan {plan}", flush=True)
    if plan in (4, 5, 6):
        s.set_angular(1)
    if plan in (0, 4, 5):
        ref = d.rhs(u0, H, dH, ubg, wl.gamma)
        s.set_gemm_plan(plan, 5, 1)
        one = s.rhs(dev(u0)).cpu().numpy()
        rnd = _pin_split(s, plan)
        got = s.rhs(dev(u0)).cpu().numpy()
        scale = max(np.max(np.abs(ref)), _term_scale(d, u0))
    elif plan in (1, 6):
        ref = d.apply_filter(u0)
        s.set_gemm_plan(plan, 5, 1)
        one = s.filter(dev(u0)).cpu().numpy()
        rnd = _pin_split(s, plan)
        got = s.filter(dev(u0)).cpu().numpy()
        scale = np.max(np.abs(ref))
    else:
        s.set_gemm_plan(plan, 5, 1)
        _, one = _step_dot(d, s, wl, u0, ubg, H, dH, plan)
        rnd = _pin_split(s, plan)
        err, got = _step_dot(d, s, wl, u0, ubg, H, dH, plan)
        print(f"  round, chunks {rnd}: step transpose dot test {err:.2e}", flush=True)
        assert err < 1e-12
        scale = np.max(np.abs(one))
        ref = one
    e_or = np.max(np.abs(got - ref)) / scale
    e_one = np.max(np.abs(got - one)) / scale
    print(f"  round, chunks {rnd}: vs oracle {e_or:.2e}, vs one launch {e_one:.2e}", flush=True)
    assert e_or < 1e-12 and e_one < 1e-13
    s.close()


@pytest.mark.parametrize("plan", [7, 8, 9, 10])
def test_split_plans_of_the_tensor_filter(plan):
    params = (2.0 / 3.0, 36.0, 8.0)
    wl, d, s, u0, ubg, H, dH = _setup(2, params)
    print(f"\n[case] forced split of GEMM plan {plan} (tensor-coupled filter)", flush=True)
    if plan in (7, 8):
        ref = d.apply_filter(u0)
        s.set_gemm_plan(plan, 5, 1)
        one = s.filter(dev(u0)).cpu().numpy()
        rnd = _pin_split(s, plan)
        got = s.filter(dev(u0)).cpu().numpy()
        scale = np.max(np.abs(ref))
    else:
        s.set_gemm_plan(plan, 5, 1)
        _, one = _step_dot(d, s, wl, u0, ubg, H, dH, plan)
        rnd = _pin_split(s, plan)
        err, got = _step_dot(d, s, wl, u0, ubg, H, dH, plan)
        print(f"  round, chunks {rnd}: step transpose dot test {err:.2e}", flush=True)
        assert err < 1e-12
        ref = one
        scale = np.max(np.abs(one))
    e_or = np.max(np.abs(got - ref)) / scale
    e_one = np.max(np.abs(got - one)) / scale
    print(f"  round, chunks {rnd}: vs oracle {e_or:.2e}, vs one launch {e_one:.2e}", flush=True)
    assert e_or < 1e-12 and e_one < 1e-13
    s.close()


def test_pinning_rejects_bad_plans():
    wl, d, s, u0, ubg, H, dH = _setup(0, None)
    for args in ((11, 5, 1, -1, 0, 0), (1, 5, 1, -1, 0, 0), (4, 5, 1, -1, 0, 0), (0, 5, 3, -1, 0, 0),
                 (0, 5, 1, 0, 9, 4), (0, 5, 1, 0, 2, -1)):
        with pytest.raises(ghmi.GHError):
            s.set_gemm_plan(*args)
    s.set_gemm_plan(0, 5, 1)
    assert s.query(6) == 5 and s.query(14) == -1
    s.close()

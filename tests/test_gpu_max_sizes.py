"""The largest shells the library accepts, against the oracle through the C
interface: L = 63 (S = 8192 points per sphere, dense angular operators of
8192 x 16384, the 64-row theta kernel of the transform method) and n_r = 256
(the point form of the radial derivative, the column kernel's registers being
sized for fewer points).

Bars.  Every FP64 evaluation of a derivative carries a rounding error of
order eps times kappa = max(|D_r| |u| + |Theta| |u| / r + |Phi| |u| / (r sin theta))
(the standard bound for a sum of products; the operators traced from the
oracle's transforms).  kappa grows with the operator norms, like L^2 and
n_r^2: at L = 63 it is about 1e3 times the term scale, and the two sides
differ by 2.6e-12 of the term scale, above the 1e-12 the smaller tests meet.
So the RHS is compared at 1e-14 kappa (about 45 ulps of it), five steps at
n_r = 256 at the sum of those errors times dt plus the filter's roundoff, and
the filter, a product with entries of size 1, at 1e-12 of the state."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi  # noqa: E402
from parity_util import rounding_scale, rounding_scale_by_shifts  # noqa: E402
from test_gpu_parity import Case, _wl, dev  # noqa: E402

pytestmark = pytest.mark.gpu

MILD = (0.5, 0.1, 2.0)


def _kappa(c, u):
    return max(rounding_scale(c.d, j, b) for j, b in enumerate(c.d.split(u, 50)))


def _rhs_error(c, label, ref, scale):
    got = c.s.rhs(dev(c.u0)).cpu().numpy()
    diff = np.max(np.abs(got - ref))
    print(f"  {label}: rhs max diff {diff:.3e}, / scale {scale:.3e} = {diff / scale:.3e}", flush=True)
    return diff / scale


@pytest.fixture(scope="module")
def deg63():
    """One shell of the largest degree: the library context (host operators of
    8192 x 16384 built and tuned) and the oracle domain; the oracle's RHS and
    rounding scale are added by the first test that needs them."""
    import time
    t0 = time.perf_counter()
    wl = _wl("L63", [(0, 3, 63, 1.8, 2.2)], [(1.0, 0.3, (0.2, 0.3, 0.4))], dt=[1e-4], filt=configs.FILTER_DEFAULT)
    c = Case(wl, pert_amp=1e-3, seed=21)
    print(f"  L = 63 context, oracle domain and inputs ready in {time.perf_counter() - t0:.1f} s", flush=True)
    return {"c": c}


def _oracle63(st, what):
    """The oracle's RHS, rounding scale or filtered state of the L = 63 case,
    each computed once (about 10 to 20 s of host time each)."""
    c = st["c"]
    if what not in st:
        if what == "ref":
            st[what] = c.oracle_rhs(c.u0)
        elif what == "kappa":
            st[what] = rounding_scale_by_shifts(c.d, 0, c.d.split(c.u0, 50)[0])
        else:
            st[what] = c.d.apply_filter(c.u0)
    return st[what]


def test_largest_degree_context(deg63):
    c = deg63["c"]
    assert c.s.P == 3 * 8192 and c.s.query(8) == 0


@pytest.mark.parametrize("what", ["ref", "kappa", "fref"])
def test_largest_degree_oracle(deg63, what):
    v = np.asarray(_oracle63(deg63, what))
    assert np.all(np.isfinite(v)) and np.max(np.abs(v)) > 0


def test_largest_degree_dense(deg63):
    c = deg63["c"]
    ref, kappa, fref = (_oracle63(deg63, w) for w in ("ref", "kappa", "fref"))
    assert _rhs_error(c, "L = 63 dense (scale kappa)", ref, kappa) < 1e-14
    got = c.s.filter(dev(c.u0)).cpu().numpy()
    ef = np.max(np.abs(got - fref)) / np.max(np.abs(fref))
    print(f"  L = 63 exponential filter: rel err {ef:.3e}", flush=True)
    assert ef < 1e-12


def test_largest_degree_by_transforms(deg63):
    c = deg63["c"]
    ref, kappa, fref = (_oracle63(deg63, w) for w in ("ref", "kappa", "fref"))
    c.s.set_angular(1)
    assert c.s.query(9) == 1 and c.s.query(10) == 1
    assert _rhs_error(c, "L = 63 by transforms (scale kappa)", ref, kappa) < 1e-14
    got = c.s.filter(dev(c.u0)).cpu().numpy()
    ef = np.max(np.abs(got - fref)) / np.max(np.abs(fref))
    print(f"  L = 63 filter by transforms: rel err {ef:.3e}", flush=True)
    assert ef < 1e-12
    c.s.set_angular(0)


def test_most_radial_points():
    rmin = configs.min_radial_spacing(256, 1.8, 2.2)
    wl = _wl("nr256", [(0, 256, 3, 1.8, 2.2)], [(1.0, 0.3, (0.2, 0.3, 0.4))], dt=[0.25 * rmin], filt=MILD)
    c = Case(wl, pert_amp=1e-3, seed=22)
    kappa = _kappa(c, c.u0)
    assert _rhs_error(c, "n_r = 256 (scale kappa)", c.oracle_rhs(c.u0), kappa) < 1e-14
    u = dev(c.u0)
    c.s.step(u, 5)
    ref = c.u0.copy()
    for _ in range(5):
        ref = c.d.rk3_step(ref, c.H, c.dH, c.ubg, c.wl.gamma, c.wl.dt)
    got = u.cpu().numpy()
    # each stage adds dt times an RHS error below 1e-14 kappa, and the filter
    # acts on O(1) data with roundoff below 1e-14 of the state
    bound = 5 * (wl.dt[0] * 1e-14 * kappa + 1e-14 * np.max(np.abs(ref)))
    diff = np.max(np.abs(got - ref))
    print(f"  5 steps: max diff {diff:.3e}, bound {bound:.3e}, change {np.max(np.abs(ref - c.u0)):.3e}",
          flush=True)
    assert diff < bound

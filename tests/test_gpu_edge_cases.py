"""Edge cases of the path against the oracle, through the C interface.

* the smallest shells the library accepts (n_r = 3, L = 1: S = 8, a 150 x 16
  x 8 GEMM far below every tile) next to a large-L instance, with a mild
  filter (the default one would remove every l = 1 degree of the metric at
  L = 1, and the evolution then loses its Lorentzian metric after one step,
  in the oracle as on the GPU);
* the exact Kerr-Schild state with no perturbation (the RHS is pure
  truncation error, a near-cancellation of large terms);
* zero steps leave the state bitwise unchanged; a negative count, a null or
  aliased pointer and an unknown kernel kind are errors;
* the transform method and the tensor-coupled filter at L = 1.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import domain  # noqa: E402
from paper_1804_09101_amd import configs, ghmi  # noqa: E402
from test_gpu_parity import Case, _wl, dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _check_rhs(c, u0, label):
    got = c.s.rhs(dev(u0)).cpu().numpy()
    ref = c.oracle_rhs(u0)
    scale = max(np.max(np.abs(ref)), c.term_scale(u0))
    err = np.max(np.abs(got - ref)) / scale
    print(f"  {label}: rhs rel err {err:.3e}", flush=True)
    assert err < 1e-12


def test_smallest_shells_next_to_a_large_instance():
    shells = [(0, 3, 1, 1.8, 2.2), (0, 3, 1, 2.2, 2.9), (1, 5, 11, 1.7, 3.0)]
    holes = [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0.3, -0.2, 0.9))]
    wl = _wl("smallest", shells, holes, filt=(0.5, 0.1, 2.0))
    c = Case(wl, pert_amp=1e-3, seed=11)
    _check_rhs(c, c.u0, "n_r = 3, L = 1 next to L = 11")
    u = dev(c.u0)
    c.s.step(u, 10)
    ref = c.u0.copy()
    for _ in range(10):
        ref = c.d.rk3_step(ref, c.H, c.dH, c.ubg, c.wl.gamma, c.wl.dt)
    err = np.max(np.abs(u.cpu().numpy() - ref)) / np.max(np.abs(ref - c.u0))
    print(f"  10 filtered steps: err/change {err:.3e}", flush=True)
    assert err < 1e-10
    c.s.set_angular(1)
    _check_rhs(c, c.u0, "L = 1 by transforms")


def test_exact_kerr_schild_state():
    wl = _wl("exact_ks", [(0, 9, 7, 1.8, 3.0), (0, 9, 7, 3.0, 5.0)], [(1.0, 0.6, (0.2, 0.3, 0.4))])
    c = Case(wl, pert_amp=0.0)
    _check_rhs(c, c.u0, "exact Kerr-Schild")


def test_tensor_filter_at_L1():
    shells = [(0, 3, 1, 1.8, 2.2), (0, 4, 1, 2.2, 2.9)]
    wl = _wl("tf_L1", shells, [(1.0, 0.0, (0, 0, 1))])
    params = (0.0, 3.0, 2.0)
    d = domain.Domain([domain.Shell(*s) for s in shells], filter_params=params, filter_kind=2)
    u0, ubg, H, dH = wl.initial_data(d.xyz(), d.offsets)
    u = u0 + 1e-3 * np.random.default_rng(3).standard_normal(u0.shape)
    s = ghmi.GHSolver(shells, 1, params, filter_kind=2)
    got = s.filter(dev(u)).cpu().numpy()
    ref = d.apply_filter(u)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"  tensor filter at L = 1: rel err {err:.3e}", flush=True)
    assert err < 1e-12


def test_zero_steps_and_argument_errors():
    c = Case(configs.single_shell(), pert_amp=1e-3, seed=2)
    u = dev(c.u0)
    before = u.clone()
    c.s.step(u, 0)
    torch.cuda.synchronize()
    assert torch.equal(u, before)
    with pytest.raises(ghmi.GHError) as ei:
        c.s._check(c.s.lib.gh_step(c.s.h, ghmi.ctypes.c_void_p(u.data_ptr()), -1))
    assert ei.value.code == -1
    with pytest.raises(ghmi.GHError) as ei:
        c.s._check(c.s.lib.gh_rhs(c.s.h, None, ghmi.ctypes.c_void_p(u.data_ptr())))
    assert ei.value.code == -1
    with pytest.raises(ghmi.GHError) as ei:
        c.s._check(c.s.lib.gh_rhs(c.s.h, ghmi.ctypes.c_void_p(u.data_ptr()), ghmi.ctypes.c_void_p(u.data_ptr())))
    assert ei.value.code == -1
    n = ghmi.ctypes.c_longlong()
    ms = ghmi.ctypes.c_double()
    with pytest.raises(ghmi.GHError) as ei:
        c.s._check(c.s.lib.gh_kernel_stats(c.s.h, len(ghmi.KERNEL_KINDS), ghmi.ctypes.byref(n), ghmi.ctypes.byref(ms)))
    assert ei.value.code == -1

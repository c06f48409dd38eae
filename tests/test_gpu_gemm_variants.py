"""Every kernel variant of the grouped GEMM, in every tile order, pinned in
turn (gh_set_gemm_variant) for the derivative and the filter GEMM, on a
mixed-L domain whose sizes are ragged for every tile: K = S = 72 (L = 5, not a
multiple of 16 or 32), 128 and 288; row counts 50 n_r not multiples of the tile
heights.  The RHS must match the oracle to 1e-12 of the term scale and a
filtered step the autotuned one to 1e-13 of the state."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_1804_09101_amd import configs, ghmi  # noqa: E402
from test_gpu_parity import Case, _wl, dev  # noqa: E402

pytestmark = pytest.mark.gpu


def test_every_variant_and_order():
    shells = [(0, 7, 5, 1.8, 2.7), (0, 9, 5, 2.7, 4.0), (1, 5, 7, 1.7, 2.9), (2, 6, 11, 1.6, 3.1)]
    holes = [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0.3, -0.2, 0.9)), (0.9, 0.2, (0.1, 0.1, 1.0))]
    wl = _wl("variants", shells, holes, filt=configs.FILTER_DEFAULT)
    c = Case(wl, pert_amp=1e-3, seed=9)
    u = dev(c.u0)
    ref = c.oracle_rhs(c.u0)
    scale = max(np.max(np.abs(ref)), c.term_scale(c.u0))
    tuned = u.clone()
    c.s.step(tuned, 1)
    worst_rhs = worst_step = 0.0
    for shape in range(ghmi.NUM_GEMM_VARIANTS):
        for order in (0, 1, 2):
            c.s.set_gemm_variant(0, shape, order)
            c.s.set_gemm_variant(1, shape, order)
            assert c.s.query(6) == shape and c.s.query(7) == shape and c.s.query(4) == order
            got = c.s.rhs(u).cpu().numpy()
            e = np.max(np.abs(got - ref)) / scale
            v = u.clone()
            c.s.step(v, 1)
            es = float((v - tuned).abs().max() / tuned.abs().max())
            print(f"  variant {shape} order {order}: rhs {e:.2e}, filtered step vs tuned {es:.2e}", flush=True)
            worst_rhs, worst_step = max(worst_rhs, e), max(worst_step, es)
            assert e < 1e-12 and es < 1e-13
    for bad in ((2, 0, 0), (0, ghmi.NUM_GEMM_VARIANTS, 0), (0, 0, 3), (0, -1, 0)):
        with pytest.raises(ghmi.GHError) as ei:
            c.s.set_gemm_variant(*bad)
        assert ei.value.code == -1


def test_misaligned_state_runs_on_the_staged_twin():
    """The direct-to-LDS variants (13-16) move A with 16-byte loads; a state
    whose base is only 8-byte aligned (a view one double into a buffer) runs on
    the register-staged twin of the same tile, which accumulates in the same
    order: bitwise the same RHS, and the oracle's to 1e-12."""
    shells = [(0, 7, 7, 1.8, 2.7), (0, 9, 7, 2.7, 4.0), (1, 6, 11, 1.6, 3.1)]
    holes = [(1.0, 0.0, (0, 0, 1)), (1.0, 0.5, (0.3, -0.2, 0.9))]
    c = Case(_wl("misaligned", shells, holes), pert_amp=1e-3, seed=5)
    u = dev(c.u0)
    buf = torch.empty(u.numel() + 1, dtype=torch.float64, device=u.device)
    um = buf[1:]
    um.copy_(u)
    assert u.data_ptr() % 16 == 0 and um.data_ptr() % 16 == 8
    ref = c.oracle_rhs(c.u0)
    scale = max(np.max(np.abs(ref)), c.term_scale(c.u0))
    for shape in (13, 14, 15, 16, 17):
        c.s.set_gemm_variant(0, shape, 1)
        a = c.s.rhs(u)
        b = c.s.rhs(um)
        e = float(np.max(np.abs(b.cpu().numpy() - ref)) / scale)
        print(f"  variant {shape}: misaligned vs aligned {'bitwise' if torch.equal(a, b) else 'DIFFERENT'}, "
              f"vs oracle {e:.2e}", flush=True)
        assert torch.equal(a, b) and e < 1e-12


def test_split_plan_matches_one_launch():
    """pulse_8shell's derivative GEMM has 1 056 tiles of 128 x 64, 4.125 per
    CU of the MI355X: the tuner may split it into whole rounds plus a tail over
    K chunks.  Whatever it keeps, the RHS matches the oracle, and the RHS and a
    filtered step match the same variants pinned as one launch up to the
    rounding of the reordered K sums (1e-13 of the term scale and of the
    state); two runs of the split plan are bitwise equal."""
    wl = configs.pulse_8shell()
    c = Case(wl)
    u = dev(c.u0)
    tuned_rhs = c.s.rhs(u)
    assert torch.equal(c.s.rhs(u), tuned_rhs)
    tuned_step = u.clone()
    c.s.step(tuned_step, 1)
    print(f"  tuned: derivative variant {c.s.query(6)} tail {c.s.query(14)} over {c.s.query(16)} K chunks, "
          f"filter variant {c.s.query(7)} tail {c.s.query(15)}", flush=True)
    ref = c.oracle_rhs(c.u0)
    scale = max(np.max(np.abs(ref)), c.term_scale(c.u0))
    err = np.max(np.abs(tuned_rhs.cpu().numpy() - ref)) / scale
    assert err < 1e-12
    c.s.set_gemm_variant(0, c.s.query(6), c.s.query(4))
    c.s.set_gemm_variant(1, c.s.query(7), c.s.query(5))
    assert c.s.query(14) == -1 and c.s.query(15) == -1 and c.s.query(16) == 0
    one = u.clone()
    c.s.step(one, 1)
    d_rhs = float((c.s.rhs(u) - tuned_rhs).abs().max()) / scale
    d_step = float((one - tuned_step).abs().max() / one.abs().max())
    print(f"  split vs one launch: rhs {d_rhs:.2e} of the term scale, step {d_step:.2e} of the state", flush=True)
    assert d_rhs < 1e-13 and d_step < 1e-13

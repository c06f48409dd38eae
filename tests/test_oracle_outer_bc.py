"""Pins of the oracle's constraint-preserving outer boundary treatment
(gh.outer_constraint_preserving; the paper's ApplyBCs case (ii), Conclusions).

The condition is defined by what it does to the characteristic fields, so
the pins check exactly that, at random states and normals:
  * outgoing fields are untouched;
  * the incoming u^psi and u^0 no longer depend on normal derivatives: adding
    s_k w to every Cartesian derivative d_k u (any w) changes the raw d_t u,
    but not the treated incoming fields (a wrong sign, index or projector in
    the constraint terms leaves a normal-derivative dependence);
  * incoming u^- is frozen;
  * on an exact solution with exact derivatives (constraints zero) the
    treatment changes nothing but u^-;
  * on a small evolution whose pulse leaves through the outer boundary, the
    constraint norm decays with the treatment and grows with Dirichlet.
"""

import numpy as np
import pytest

from oracle import domain, gh, grid
from oracle import kerr_schild as ks
from paper_1804_09101_amd import configs, inputs


def _state(seed, npts=9):
    xyz = grid.ShellGrid(3, 2, 5.0, 6.0).xyz()[:, :npts]
    ex = ks.exact_fields(xyz, M=1.0, chi=0.6, axis=(0.2, -0.1, 1.0))
    rng = np.random.default_rng(seed)
    u = ex["u"] + 1e-2 * rng.standard_normal(ex["u"].shape)
    du = ex["du"] + 1e-2 * rng.standard_normal(ex["du"].shape)
    H = ex["H"] + 1e-3 * rng.standard_normal(ex["H"].shape)
    dH = ex["dH"].reshape(4, 4, -1)
    n = xyz / np.sqrt(np.sum(xyz * xyz, axis=0))       # outward radial normal
    return u, du, H, dH, n


def _treat(u, du, H, dH, n, gam):
    psi, _, _ = gh.unpack_fields(u)
    geo = gh.Geometry(psi)
    s_lo, s_up = gh.unit_normal(geo, n)
    raw = gh.rhs_pointwise(u, du, H, dH, *gam)
    out = gh.outer_constraint_preserving(raw, u, du, s_lo, s_up, geo, gam[1], gam[2])
    return raw, out, geo, s_lo, s_up


@pytest.mark.parametrize("gam", [(1.0, -1.0, 1.0), (0.4, 0.5, 1.3), (1.0, -0.3, 0.0)])
def test_outgoing_untouched_incoming_free_of_normal_derivatives(gam):
    u, du, H, dH, n = _state(1)
    raw, out, geo, s_lo, s_up = _treat(u, du, H, dH, n, gam)
    v_psi, v_0, v_p, v_m = gh.char_speeds(geo, s_lo, gam[1])
    assert np.all(v_0 < 0) and np.all(v_m < 0) and np.all(v_p > 0)   # outward shift at r ~ 5
    f_raw = gh.char_fields(raw, s_lo, s_up, gam[2])
    f_out = gh.char_fields(out, s_lo, s_up, gam[2])
    assert np.max(np.abs(f_out[2] - f_raw[2])) < 1e-15 * np.max(np.abs(f_raw[2]))   # u^+ untouched
    assert np.max(np.abs(f_out[3])) < 1e-15 * np.max(np.abs(f_raw[3]))                # u^- frozen
    # normal derivatives changed by s_k w
    w = np.random.default_rng(2).standard_normal((50, u.shape[1]))
    du2 = du + s_lo[:, None, :] * w[None]
    raw2, out2, _, _, _ = _treat(u, du2, H, dH, n, gam)
    f_raw2 = gh.char_fields(raw2, s_lo, s_up, gam[2])
    f_out2 = gh.char_fields(out2, s_lo, s_up, gam[2])
    assert np.max(np.abs(f_raw2[1] - f_raw[1])) > 1e-3                 # the raw u^0 does depend on them
    assert np.max(np.abs(f_out2[1] - f_out[1])) < 1e-13                # the treated u^0 does not
    incoming_psi = v_psi < 0
    if np.any(incoming_psi):
        assert np.max(np.abs(f_raw2[0] - f_raw[0])) > 1e-3
        assert np.max(np.abs((f_out2[0] - f_out[0])[:, incoming_psi])) < 1e-13
    else:
        # gamma1 = -1: u^psi has speed zero and is left as it is
        assert np.max(np.abs(f_out[0] - f_raw[0])) < 1e-15
    assert np.max(np.abs(f_out2[2] - f_raw2[2])) < 1e-14                # u^+ still the raw one


def test_exact_solution_is_left_alone_except_incoming_u_minus():
    """A boosted hole with exact derivatives: every constraint vanishes, so the
    treated u^psi and u^0 equal the exact time derivatives' projections."""
    xyz = grid.ShellGrid(3, 2, 5.0, 6.0).xyz()[:, :12]
    ex = ks.exact_fields(xyz, M=1.0, chi=0.4, axis=(0.1, 0.5, 0.3), boost=(0.2, -0.1, 0.15))
    gam = (0.7, 0.4, 1.1)
    n = xyz / np.sqrt(np.sum(xyz * xyz, axis=0))
    raw, out, geo, s_lo, s_up = _treat(ex["u"], ex["du"], ex["H"], ex["dH"].reshape(4, 4, -1), n, gam)
    assert np.max(np.abs(raw - ex["dtu"])) < 1e-13
    f_ex = gh.char_fields(ex["dtu"], s_lo, s_up, gam[2])
    f_out = gh.char_fields(out, s_lo, s_up, gam[2])
    for j in (0, 1, 2):
        assert np.max(np.abs(f_out[j] - f_ex[j])) < 1e-13
    assert np.max(np.abs(f_ex[3])) > 1e-3 and np.max(np.abs(f_out[3])) < 1e-15 * np.max(np.abs(f_ex[3]))


def test_constraint_norm_decays_with_the_treatment_and_grows_with_dirichlet():
    shells = [(0, 9, 5, 1.8, 3.5), (0, 9, 5, 3.5, 6.0)]
    wl = configs.Workload("cpbc", shells, [(1.0, 0.0, (0, 0, 1))], [(1.0, -1.0, 1.0)], [0.0125],
                          configs.FILTER_DEFAULT, 160, None)
    norms = {}
    for bc in ("dirichlet", "constraint_preserving"):
        d = domain.Domain([domain.Shell(*s) for s in shells], filter_params=configs.FILTER_DEFAULT, outer_bc=bc)
        u0, ubg, H, dH = wl.initial_data(d.xyz(), d.offsets)
        u = u0 + d.to_layout(inputs.gaussian_pulse_Pi(d.xyz(), 1e-3, 5.0, 0.5, 0))
        n0 = d.constraint_norm(u, H)[0]
        for _ in range(160):
            u = d.rk3_step(u, H, dH, ubg, wl.gamma, wl.dt)
        norms[bc] = (n0, d.constraint_norm(u, H)[0])
    (n0, nd), (_, nc) = norms["dirichlet"], norms["constraint_preserving"]
    assert nc < 0.5 * n0 and nd > 1.5 * n0 and nd > 3.0 * nc
